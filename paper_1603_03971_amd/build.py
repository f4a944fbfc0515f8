"""Build librtm.so (HIP, gfx950) in-tree with hipcc, and the stand-alone bandwidth probe.

Flags: FP contraction off (the kernels spell out every FMA, so halo and interior agree bitwise),
packed-FP32 instructions off, fast hardware float atomics for injection.  The two sources compile
in parallel to objects under _build/, which are then linked into the shared library.  The probe
(csrc/stream_probe.hip, a program of its own that the library does not use) is built beside it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "rtm.hip"), os.path.join(HERE, "csrc", "cnn.hip")]
LIB = os.path.join(HERE, "librtm.so")
PROBE_SRC = os.path.join(HERE, "csrc", "stream_probe.hip")
PROBE = os.path.join(HERE, "stream_probe")
OBJDIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("RTM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-ffp-contract=off", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(os.path.basename(src))[0] + ".o")
        cmd = ["hipcc", *FLAGS, *extra, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    probe_cmd = ["hipcc", "-O3", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
                 "-packed-fp32-ops", "-o", PROBE + ".tmp", PROBE_SRC]
    procs.append((probe_cmd, subprocess.Popen(probe_cmd)))
    for cmd, p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    os.replace(PROBE + ".tmp", PROBE)
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs, "-ldl"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
