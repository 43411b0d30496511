"""Compile the gfx950 C-ABI library libwave.so in-tree with hipcc.

The step kernels of each space order are a translation unit of their own
(csrc/wave_o<order>.hip), so the units compile in parallel (at most MAX_JOBS
at once, default: the CPU count).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libwave.so")
ORDERS = (2, 4, 6, 8, 10, 12, 14, 16)
SOURCES = ["wave_host.cpp", "wave_kernels.hip"] + [f"wave_o{o}.hip" for o in ORDERS]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions; arithmetic exactly as written (explicit fmaf only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-result", "-Wno-c++20-extensions",
]


def build(verbose: bool = False, out_dir: str = OUT, defines=(), jobs: int = 0, orders=ORDERS,
          extra_flags=()) -> str:
    """Compile libwave.so into ``out_dir``.  ``defines`` and ``orders`` serve
    experimental builds (extra ``-D`` knobs; a single space order, which then
    also restricts the order dispatch)."""
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, "libwave.so")
    jobs = jobs or int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 4
    orders = tuple(orders)
    if orders != ORDERS:
        if len(orders) != 1:
            raise ValueError("an experimental build holds all orders or exactly one")
        defines = tuple(defines) + (f"WAVE_ONLY_ORDER={orders[0]}",)
    pending = ["wave_host.cpp", "wave_kernels.hip"] + [f"wave_o{o}.hip" for o in orders]
    running = []
    objs = []
    failed = []
    while pending or running:
        while pending and len(running) < jobs:
            src = pending.pop(0)
            obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
            cmd = [HIPCC, *FLAGS, *extra_flags, *[f"-D{d}" for d in defines], "-c",
                   os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                  stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        src, proc = running.pop(0)
        out, _ = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(out)
            failed.append(src)
        elif verbose:
            warn = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
            if warn:
                print("\n".join(warn), flush=True)
    if failed:
        raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
