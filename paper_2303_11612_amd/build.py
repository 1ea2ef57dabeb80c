"""Build the HIP library in-tree for gfx950.

``python -m paper_2303_11612_amd.build`` (or ``build()``) compiles the
translation units under ``csrc/`` (in parallel) and links them into
``libtucker_rand.so`` next to this file.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# translation units, compiled in parallel and linked into one library: the
# host driver, the factor kernel instances, the low-precision power steps and
# the batched driver
SOURCES = [
    # one unit per factor kernel instance (FactorVariant 0 .. 15), the slowest
    ("tr_factor_inst.hip", (f"-DTR_FACTOR_INST={k}",)) for k in range(17)] + [
    ("tr_lowp_launch.hip", ()), ("tucker_rand.hip", ()), ("tr_factor_launch.hip", ()),
    ("tr_pw_fused.hip", ()), ("tr_batch.hip", ())]
SRC = os.path.join(CSRC, "tucker_rand.hip")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtucker_rand.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False, extra_flags=()) -> str:
    import tempfile
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="tucker_rand_build_") as tmpdir:
        objs, cmds = [], []
        for k, (src, defs) in enumerate(SOURCES):
            obj = os.path.join(tmpdir, f"{k:02d}_" + os.path.splitext(src)[0] + ".o")
            cmds.append((src, [cc, *HIPCC_FLAGS, *defs, *extra_flags, "-I", INCLUDE, "-I", CSRC,
                               "-c", os.path.join(CSRC, src), "-o", obj]))
            objs.append(obj)
        # the factor instances dominate; run them first, at most one per core
        jobs = max(1, min(len(cmds), os.cpu_count() or 1))
        failed, running, queue = [], [], list(reversed(cmds))
        while queue or running:
            while queue and len(running) < jobs:
                src, cmd = queue.pop()
                if verbose:
                    print(" ".join(cmd), flush=True)
                running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                      stderr=subprocess.STDOUT, text=True)))
            src, pr = running.pop(0)
            out, _ = pr.communicate()
            if pr.returncode != 0:
                failed.append((src, out))
            elif verbose and out.strip():
                sys.stderr.write(out)
        if failed:
            for src, out in failed:
                sys.stderr.write(f"--- {src}\n{out}")
            raise RuntimeError(f"hipcc failed for {', '.join(s for s, _ in failed)}")
        tmp = LIB + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"link failed with exit code {res.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
