"""Build the host-sanitizer driver: a copy of libhfx.so whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer (device code as in the main
build, whose objects are reused), and hostsan_driver linked against it with
the sanitizer runtime inside the executable.  Output: tests/hostsan/_build/."""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
MAIN = os.path.join(ROOT, "paper_2009_03559_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build():
    os.makedirs(OUT, exist_ok=True)
    for d in ("gen", "obj"):
        src, dst = os.path.join(MAIN, d), os.path.join(OUT, d)
        if os.path.isdir(src) and not os.path.isdir(dst):
            shutil.copytree(src, dst)
    env = dict(os.environ, HFX_BUILD_DIR=OUT, HFX_HOST_SANITIZE="1")
    subprocess.check_call([sys.executable, os.path.join(ROOT, "paper_2009_03559_amd", "build.py"), "--changed"],
                          env=env)
    exe = os.path.join(OUT, "hostsan_driver")
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17"] + SAN +
                          ["-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "hostsan_driver.cpp"),
                           "-o", exe, "-L" + OUT, "-lhfx", "-Wl,-rpath," + OUT])
    return exe


if __name__ == "__main__":
    print(build())
