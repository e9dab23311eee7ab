"""Build the test helper librocrand_probe.so (host-only use of rocRAND's
Philox4x32-10 engine, an external reference for the Philox pins)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librocrand_probe.so")


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.check_call(
        ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-fPIC", "-shared", "-x", "hip",
         os.path.join(HERE, "rocrand_probe.cpp"), "-o", tmp],
        stderr=subprocess.DEVNULL)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
