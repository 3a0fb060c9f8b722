"""Builds the plain C client of librtm (rtm_c_demo) next to its source: gcc,
the public header and the HIP runtime only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))


def build() -> str:
    out = os.path.join(HERE, "rtm_c_demo")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
           os.path.join(HERE, "rtm_c_demo.c"),
           "-L" + os.path.join(ROOT, "paper_2201_06914_amd"), "-lrtm",
           "-L/opt/rocm/lib", "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_2201_06914_amd", "-Wl,-rpath,/opt/rocm/lib",
           "-o", out]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build())
