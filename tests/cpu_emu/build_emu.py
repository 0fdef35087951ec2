"""Build the library's kernel sources as a CPU program (see hip/hip_runtime.h here)."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2207_04649_amd", "csrc")


def build(out_dir: str, asan: bool = False, defines: tuple = ()) -> str:
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
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(tmp, exe)
    return exe
