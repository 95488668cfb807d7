"""Build libnegf_hostsim.so: the library's host orchestration (csrc/api.hip)
linked with the CPU test double of its kernels (hostsim.cpp).  CPU tests only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2602_03438_amd", "csrc")
LIB = os.path.join(HERE, "libnegf_hostsim.so")


LIB_SANITIZED = os.path.join(HERE, "libnegf_hostsim_sanitized.so")
# host code only: AddressSanitizer and UndefinedBehaviorSanitizer (every finding fatal)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """The shared AddressSanitizer runtime of the compiler that builds the sanitized library (a
    process that loads the library must preload it)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    r = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], check=True, capture_output=True,
                       text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path):
        r = subprocess.run([hipcc, "-print-resource-dir"], check=True, capture_output=True, text=True)
        path = os.path.join(r.stdout.strip(), "lib", "linux", "libclang_rt.asan-x86_64.so")
    return path


def build(sanitize: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = os.path.join(ROOT, "_build", "hostsim_sanitized" if sanitize else "hostsim")
    os.makedirs(out, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-Wno-unused-result"] + (SANITIZE if sanitize else [])
    objs = []
    for src in (os.path.join(CSRC, "api.hip"), os.path.join(CSRC, "serinv.hip"), os.path.join(HERE, "hostsim.cpp")):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        subprocess.run([hipcc, *flags, "-x", "hip", "-c", src, "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    lib = LIB_SANITIZED if sanitize else LIB
    link = ["-shared-libasan", *SANITIZE] if sanitize else []
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *link, "-o", lib, *objs], check=True,
                   capture_output=True)
    return lib


if __name__ == "__main__":
    import sys
    print(build(sanitize="--sanitize" in sys.argv))
