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


LIB_TSAN = os.path.join(HERE, "libnegf_hostsim_tsan.so")
# host code only: ThreadSanitizer
SANITIZE_THREAD = ["-Xarch_host", "-fsanitize=thread", "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime(name: str = "asan") -> str:
    """The shared sanitizer runtime (``asan`` or ``tsan``) of the compiler that builds the
    sanitized library (a process that loads the library must preload it)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = f"libclang_rt.{name}-x86_64.so"
    r = subprocess.run([hipcc, f"-print-file-name={lib}"], check=True, capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path):
        r = subprocess.run([hipcc, "-print-resource-dir"], check=True, capture_output=True, text=True)
        path = os.path.join(r.stdout.strip(), "lib", "linux", lib)
    return path


def asan_runtime() -> str:
    return runtime("asan")


def build(sanitize=False) -> str:
    """sanitize: False, True (AddressSanitizer + UndefinedBehaviorSanitizer) or "thread"."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tsan = sanitize == "thread"
    out = os.path.join(ROOT, "_build", "hostsim_tsan" if tsan else "hostsim_sanitized" if sanitize else "hostsim")
    os.makedirs(out, exist_ok=True)
    san = SANITIZE_THREAD if tsan else SANITIZE if sanitize else []
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-Wno-unused-result"] + san
    objs = []
    for src in (os.path.join(CSRC, "api.hip"), os.path.join(CSRC, "serinv.hip"), os.path.join(HERE, "hostsim.cpp")):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        subprocess.run([hipcc, *flags, "-x", "hip", "-c", src, "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    lib = LIB_TSAN if tsan else LIB_SANITIZED if sanitize else LIB
    link = SANITIZE_THREAD if tsan else ["-shared-libasan", *SANITIZE] if sanitize else []
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *link, "-o", lib, *objs], check=True,
                   capture_output=True)
    return lib


if __name__ == "__main__":
    import sys
    print(build(sanitize="thread" if "--tsan" in sys.argv else "--sanitize" in sys.argv))
