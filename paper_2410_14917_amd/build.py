"""Build libkrylov_phi.so in-tree with hipcc for gfx950, and the C-ABI test
client (tests/c_abi_client: host C++ against the HIP runtime and the library,
no Python)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "krylov_phi.hip")
OUT = os.path.join(HERE, "libkrylov_phi.so")
TIMELINE_OUT = os.path.join(HERE, "libkrylov_phi_timeline.so")
CLIENT_SRC = os.path.join(ROOT, "tests", "c_abi_client.cpp")
CLIENT = os.path.join(ROOT, "tests", "c_abi_client")
RUNNER_SRC = os.path.join(HERE, "kp_run.cpp")
RUNNER = os.path.join(HERE, "kp_run")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    cmd = [hipcc, *FLAGS, SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, OUT)
    build_timeline(verbose)
    build_client(verbose)
    build_runner(verbose)
    return OUT


def build_timeline(verbose: bool = False) -> str:
    """The same library with the device timeline compiled in (KP_TIMELINE:
    kp_set_timeline records per-phase clock stamps), for profiling only."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = TIMELINE_OUT + ".tmp"
    cmd = [hipcc, *FLAGS, "-DKP_TIMELINE", SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc (timeline build) failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, TIMELINE_OUT)
    return TIMELINE_OUT


def build_runner(verbose: bool = False) -> str:
    """The native runner (kp_run.cpp: the C ABI and the system HIP runtime,
    for profiling a process that maps one runtime), next to the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = RUNNER + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), RUNNER_SRC, "-o", tmp, "-L" + HERE,
           "-lkrylov_phi", "-Wl,-rpath,$ORIGIN"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("building kp_run failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, RUNNER)
    return RUNNER


def build_client(verbose: bool = False) -> str:
    """Host-only program: g++ with the HIP runtime headers; it finds the
    library next to it in the tree through an $ORIGIN-relative rpath."""
    cxx = os.environ.get("CXX", "g++")
    tmp = CLIENT + ".tmp"
    cmd = [cxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROCM, "include"), CLIENT_SRC, "-o", tmp, "-L" + HERE,
           "-lkrylov_phi", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../paper_2410_14917_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("building the C-ABI client failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, CLIENT)
    return CLIENT


if __name__ == "__main__":
    print(build(verbose=True))
