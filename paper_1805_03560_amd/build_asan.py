"""Host-side sanitizer build of the library's host code (test infrastructure).

Compiles every csrc/*.hip translation unit for the host only (no device code) with
AddressSanitizer and UndefinedBehaviorSanitizer, adds the driver tests/asan/host_checks.cpp and
links the executable _build/asan/whmc_host_checks with the clang sanitizer runtimes.  Without
device code the objects name device-image symbols that no object defines; the link gets empty
stand-ins for them, so the executable registers no usable GPU code and must not launch kernels:
the driver exercises the coefficient generators and the argument checks of every entry point,
which run before any device work.  It runs on a machine without a GPU.  Used by
tests/test_host_sanitizers.py.
"""
import concurrent.futures
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build", "asan")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
       "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
INC = ["-I", os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd[:3])} ... failed:\n{r.stderr[-6000:]}")


def _compile(src):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    _run([HIPCC, "--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950"] + SAN + INC +
         ["-c", src, "-o", obj])
    return obj


def build(jobs=None):
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with concurrent.futures.ThreadPoolExecutor(jobs or min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, srcs))
    drv = os.path.join(OUT, "host_checks.o")
    sanitize = "-fsanitize=" + "address,undefined"
    _run([CLANGXX, "-O1", "-g", "-std=c++17", sanitize, "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"] + INC +
         ["-c", os.path.join(ROOT, "tests", "asan", "host_checks.cpp"), "-o", drv])
    # empty stand-ins for the device images the host-only objects refer to
    missing = set()
    for o in objs:
        out = subprocess.run(["nm", o], capture_output=True, text=True).stdout
        missing |= {ln.split()[-1] for ln in out.splitlines() if ln.strip().startswith("U __hip_fatbin_")}
    stub_c = os.path.join(OUT, "device_image_stubs.c")
    with open(stub_c, "w") as f:
        f.write("/* generated: no device code in the host-only sanitizer build */\n")
        for name in sorted(missing):
            f.write(f"const unsigned char {name}[64] = {{0}};\n")
    stub_o = os.path.join(OUT, "device_image_stubs.o")
    _run([CLANGXX, "-x", "c", "-c", stub_c, "-o", stub_o])
    exe = os.path.join(OUT, "whmc_host_checks")
    _run([CLANGXX, sanitize, "-o", exe, drv, stub_o] + objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"])
    return exe


if __name__ == "__main__":
    print(build())
