"""Builds libcoot_front_end_cases.so, the C++ front-end test cases the GPU
tests call through ctypes (host code only: g++ against include/coot.hpp and
the library)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIBDIR = os.path.join(ROOT, "paper_2308_03120_amd")
OUT = os.path.join(HERE, "libcoot_front_end_cases.so")


def build() -> str:
    tmp = OUT + f".tmp{os.getpid()}"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", "-fPIC", "-shared",
                           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
                           os.path.join(HERE, "front_end_cases.cpp"), "-o", tmp, "-L" + LIBDIR, "-lcoot_mi355x",
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,$ORIGIN/../../paper_2308_03120_amd"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
