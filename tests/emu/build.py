"""Build the CPU emulation of libara (test infrastructure).

The library's own sources (paper_1310_2274_amd/csrc/*.hip) are compiled as
host C++ against the emulated HIP runtime in this directory, with a
sanitizer, and linked with a small driver into one executable:

    python tests/emu/build.py address|thread [out]

Every GPU thread becomes a host thread (see hip/hip_runtime.h), so
AddressSanitizer checks every device and LDS access and ThreadSanitizer
reports any cross-lane LDS access that no wave_sync / __syncthreads orders.
Host compiler only: no GPU code is built here.
"""
import fcntl
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1310_2274_amd", "csrc")
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")


def build(sanitizer: str, out: str = "") -> str:
    """Compile and link the driver; safe to call from several processes at
    once (pytest-xdist workers): one build per output at a time, objects in
    a private directory, and the executable replaced in one rename."""
    assert sanitizer in ("address", "thread")
    out = out or os.path.join(HERE, f"emu_driver_{sanitizer}")
    srcs = [os.path.join(CSRC, f) for f in ("ara_api.hip", "ara_kernels.hip", "ara_surrogate.hip")]
    cmd = [CXX, "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={sanitizer}",
           "-Wno-unknown-attributes", "-Wno-ignored-attributes", "-Wno-unused-result",
           "-I", HERE, "-I", os.path.join(ROOT, "include"), "-pthread"]
    with open(out + ".lock", "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        with tempfile.TemporaryDirectory(dir=os.path.dirname(out)) as tmp:
            objs = []
            for s in srcs + [os.path.join(HERE, "emu_runtime.cpp"), os.path.join(HERE, "emu_driver.cpp")]:
                o = os.path.join(tmp, os.path.basename(s) + ".o")
                subprocess.check_call(cmd + ["-x", "c++", "-c", s, "-o", o])
                objs.append(o)
            exe = os.path.join(tmp, "driver")
            subprocess.check_call([CXX, f"-fsanitize={sanitizer}", "-pthread", "-o", exe] + objs)
            os.replace(exe, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else "address", sys.argv[2] if len(sys.argv) > 2 else ""))
