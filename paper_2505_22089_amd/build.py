"""Build libchm.so (HIP for gfx950) in-tree, beside this file.

hipcc compiles every source of csrc/ with -O3 for gfx950 only; packed fp32
instructions are disabled for device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libchm.so")
SOURCES = ["chm_host.cpp", "sched.cpp", "driver.cpp", "sao.cpp", "ransac.cpp", "sao_device.hip", "ransac_device.hip", "project.hip", "bucket.hip", "match.hip", "match_bm.hip",
           "bruteforce.hip"]
ARCH = "gfx950"


def build(verbose: bool = False, jobs: int = 6) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["hipcc", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
              "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wall", "-Wno-unused-result"]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = common + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait() if procs[0][1].poll() is None else None
            import time
            time.sleep(0.05)
    errors = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            errors.append("%s:\n%s" % (src, text))
        elif verbose and text.strip():
            print(text)
    if errors:
        raise RuntimeError("libchm build failed:\n" + "\n".join(errors))
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print("built", OUT)
