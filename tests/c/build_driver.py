"""Compile tests/c/lb_c_driver and tests/c/lb3_c_driver (plain C programs that
drive liblb.so through include/lb.h and include/lb3.h) with gcc; run as a
script or call build()."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "lb_c_driver.c")
EXE = os.path.join(HERE, "lb_c_driver")
SRC3 = os.path.join(HERE, "lb3_c_driver.c")
EXE3 = os.path.join(HERE, "lb3_c_driver")
LIBDIR = os.path.join(ROOT, "paper_2101_04847_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def command(out: str = EXE, src: str = SRC) -> list:
    return ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), src, "-o", out,
            "-L", LIBDIR, "-llb", "-Wl,-rpath,$ORIGIN/../../paper_2101_04847_amd",
            "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]


def build(out: str = EXE, src: str = SRC) -> str:
    """Needs liblb.so built first; returns the path of the program (the 2D
    driver by default)."""
    if not os.path.exists(os.path.join(LIBDIR, "liblb.so")):
        raise RuntimeError("liblb.so is not built")
    r = subprocess.run(command(out, src), capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed building " + os.path.basename(src) + ":\n" + r.stderr)
    return out


def build_all() -> list:
    return [build(EXE, SRC), build(EXE3, SRC3)]


if __name__ == "__main__":
    print(build_all() if len(sys.argv) == 1 else build(sys.argv[1]))
