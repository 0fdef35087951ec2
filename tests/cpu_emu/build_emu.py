"""Build the library's kernel sources as a CPU program (see hip/hip_runtime.h here)."""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2207_04649_amd", "csrc")


def _stamp(cmd: list) -> str:
    """A hash of the command and of every source it reads (kernels, headers, driver)."""
    h = hashlib.sha256(" ".join(cmd).encode())
    files = sorted(glob.glob(os.path.join(CSRC, "*")) + glob.glob(os.path.join(HERE, "*.cpp")) +
                   glob.glob(os.path.join(HERE, "hip", "*")) + glob.glob(os.path.join(ROOT, "include", "*.h")))
    for f in files:
        if os.path.isfile(f):
            with open(f, "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()


def build(out_dir: str, asan: bool = False, defines: tuple = ()) -> str:
    """Builds the emulator, or reuses the one built from the same sources and options."""
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "dpc_emu_asan" if asan else "dpc_emu")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    # built under a private name and renamed into place, so that test processes
    # running side by side never execute a half-written file
    tmp = f"{exe}.{os.getpid()}.tmp"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-x", "c++", "-I", HERE, "-I", os.path.join(ROOT, "include"), *srcs,
           "-x", "none", os.path.join(HERE, "driver.cpp"), "-o", tmp]
    if asan:
        cmd[1:1] = ["-fsanitize=address", "-fno-omit-frame-pointer"]
    # extra -D options of the kernel sources (space-separated), e.g. to check a
    # compile-time variant of a kernel
    cmd[1:1] = list(defines) + os.environ.get("DPC_EMU_DEFINES", "").split()
    stamp = _stamp([c for c in cmd if c != tmp])
    stamp_file = exe + ".stamp"
    if os.path.exists(exe) and os.path.exists(stamp_file) and open(stamp_file).read() == stamp:
        return exe
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(tmp, exe)
    with open(stamp_file + f".{os.getpid()}", "w") as f:
        f.write(stamp)
    os.replace(stamp_file + f".{os.getpid()}", stamp_file)
    return exe
