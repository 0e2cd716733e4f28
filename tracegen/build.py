"""Build the trace generator libraries in-tree (host: gcc, device: hipcc)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> None:
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                    os.path.join(HERE, "tg_host.c"), "-o", os.path.join(HERE, "libtracegen_host.so")],
                   check=True)
    subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Wno-unused-result", "-Wno-unused-value",
                    os.path.join(HERE, "tg_dev.hip"), "-o", os.path.join(HERE, "libtracegen_dev.so")],
                   check=True, capture_output=True)


if __name__ == "__main__":
    build()
