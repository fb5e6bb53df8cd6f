"""Build the HIP library libnvp.so for gfx950 (hipcc; one translation unit per FFT length).

Usage: python -m paper_2011_03009_amd.build [--incremental] [-j N]
"""

import argparse
import concurrent.futures as cf
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB_DIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIB_DIR, "libnvp.so")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled: plain float code only.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE] + DEVICE_FLAGS


def lengths():
    src = open(os.path.join(CSRC, "launch.hpp")).read()
    m = re.search(r"#define NVP_FOR_EACH_LENGTH\(X\)(.*?)\n\n", src, re.S)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def _deps(src, seen=None):
    """src and the local headers it includes, transitively (quoted #include lines)."""
    seen = set() if seen is None else seen
    if src in seen or not os.path.exists(src):
        return seen
    seen.add(src)
    for inc in re.findall(r'^\s*#\s*include\s+"([^"]+)"', open(src).read(), re.M):
        _deps(os.path.normpath(os.path.join(os.path.dirname(src), inc)), seen)
    return seen


def _stale(obj, srcs):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(s) > t for s in srcs)


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build step failed: %s\n%s" % (" ".join(cmd), out))
    return out


def jobs_list():
    jobs = []
    inst = os.path.join(CSRC, "inst.hip")
    for L in lengths():
        obj = os.path.join(OBJ, "inst_%d.o" % L)
        jobs.append((obj, [HIPCC] + COMMON + ["-DNVP_L=%d" % L, "-c", inst, "-o", obj], sorted(_deps(inst))))
    for name, extra in (("kspec.hip", []), ("dispatch.cpp", []), ("runtime.cpp", ["-ffp-contract=off"]),
                        ("qbox.hip", []), ("boxnet.hip", []), ("learn.cpp", []),
                        ("incident.hip", []), ("vie.hip", []), ("noalloc.hip", []), ("difference.hip", ["-ffp-contract=off"])):
        obj = os.path.join(OBJ, os.path.splitext(name)[0] + ".o")
        jobs.append((obj, [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, name), "-o", obj],
                     sorted(_deps(os.path.join(CSRC, name)))))
    return jobs


def build(incremental=False, jobs=None, verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(LIB_DIR, exist_ok=True)
    todo = [j for j in jobs_list() if not incremental or _stale(j[0], j[2])]
    n = jobs or min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=n) as ex:
        for out in ex.map(lambda j: _run(j[1]), todo):
            if verbose and out.strip():
                print(out)
    objs = [j[0] for j in jobs_list()]
    if todo or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(incremental=a.incremental, jobs=a.j, verbose=a.v))
    sys.exit(0)
