"""Build libnegf_hostsim.so: the library's host orchestration (csrc/api.hip)
linked with the CPU test double of its kernels (hostsim.cpp).  CPU tests only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2602_03438_amd", "csrc")
LIB = os.path.join(HERE, "libnegf_hostsim.so")


def build() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = os.path.join(ROOT, "_build", "hostsim")
    os.makedirs(out, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-Wno-unused-result"]
    objs = []
    for src in (os.path.join(CSRC, "api.hip"), os.path.join(CSRC, "serinv.hip"), os.path.join(HERE, "hostsim.cpp")):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        subprocess.run([hipcc, *flags, "-x", "hip", "-c", src, "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB, *objs], check=True,
                   capture_output=True)
    return LIB


if __name__ == "__main__":
    print(build())
