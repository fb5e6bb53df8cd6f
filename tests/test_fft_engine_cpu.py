"""The Stockham FFT engine's and the source kernel's index arithmetic and synchronisation, on the CPU.

tests/fft_host/harness.cpp compiles the engine header of the library
(csrc/fft_core.hpp) for the host, runs each lane of a column as a host thread
with a barrier for every LDS exchange, and compares every use the kernels make
of it (forward with a zero upper half, inverse keeping the lower half, the
fused z-pass product with the reverse-order inverse, the even-sequence FP64
passes through the real-plane exchange, the wave-local octant-row pass, and
interleaved columns) with a direct DFT in long double, for every compiled
transform length in FP64 and FP32.  The harness is built with AddressSanitizer,
so a register or LDS index outside its array fails the test, and it checks
that every output is written exactly once.
"""

import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "fft_host")
CSRC = os.path.join(ROOT, "paper_2011_03009_amd", "csrc")
BUILD = os.path.join(HERE, "_build")


def compiled_lengths():
    src = open(os.path.join(CSRC, "launch.hpp")).read()
    m = re.search(r"#define NVP_FOR_EACH_LENGTH\(X\)(.*?)\n\n", src, re.S)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def _build_and_run(L):
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "harness_%d" % L)
    srcs = [os.path.join(HERE, "harness.cpp"), os.path.join(CSRC, "fft_core.hpp"),
            os.path.join(HERE, "hip", "hip_runtime.h")]
    if not os.path.exists(exe) or any(os.path.getmtime(s) > os.path.getmtime(exe) for s in srcs):
        cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-pthread",
               "-I" + HERE, "-I" + CSRC, "-DNVP_HOST_L=%d" % L, srcs[0], "-o", exe + ".tmp"]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            return L, False, "compile failed:\n" + r.stdout[-3000:]
        os.replace(exe + ".tmp", exe)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    return L, r.returncode == 0 and r.stdout.startswith("OK"), r.stdout[-3000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_engine_every_length_on_host_threads():
    lengths = compiled_lengths()
    assert len(lengths) >= 50 and lengths[-1] == 8192
    workers = max(1, min(8, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(_build_and_run, lengths))
    bad = [(L, out) for L, ok, out in results if not ok]
    assert not bad, "\n".join("L=%d:\n%s" % b for b in bad[:4])


def test_engine_catches_a_wrong_constant(tmp_path):
    """The harness is sharp: the same engine with one radix-9 rotation constant perturbed fails."""
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    src = open(os.path.join(CSRC, "fft_core.hpp")).read()
    bad = src.replace("0.766044443118978035202392650555", "(0.766044443118978035202392650555 + 1e-7)", 1)
    assert bad != src
    (tmp_path / "fft_core.hpp").write_text(bad)
    exe = str(tmp_path / "h")
    cmd = ["g++", "-std=c++20", "-O1", "-pthread", "-I" + HERE, "-I" + str(tmp_path), "-DNVP_HOST_L=144",
           os.path.join(HERE, "harness.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    assert r.returncode != 0 and "FAIL" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_source_kernel_on_host_threads():
    """The source kernel (csrc/source.hpp) run workgroup by workgroup on host threads against the
    transfer and source product summed directly (tests/fft_host/source_harness.cpp)."""
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "source_harness")
    srcs = [os.path.join(HERE, "source_harness.cpp"), os.path.join(CSRC, "source.hpp"),
            os.path.join(CSRC, "field_dev.hpp"), os.path.join(CSRC, "common.hpp"),
            os.path.join(CSRC, "fft_core.hpp"), os.path.join(HERE, "hip", "hip_runtime.h")]
    if not os.path.exists(exe) or any(os.path.getmtime(s) > os.path.getmtime(exe) for s in srcs):
        cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-pthread",
               "-I" + HERE, "-I" + CSRC, srcs[0], "-o", exe + ".tmp"]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, "compile failed:\n" + r.stdout[-3000:]
        os.replace(exe + ".tmp", exe)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout[-3000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_kernel_tabulation_tasks_cover_every_row_once():
    """The tasks of the kernel-tabulation pass (csrc/kz_tasks.hpp) on octant shapes of the paper's
    workloads and small edge cases: every row written once, indices in the octant, mirror pairs
    inside the square of nonzero rows (tests/fft_host/kz_tasks_check.cpp)."""
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "kz_tasks_check")
    srcs = [os.path.join(HERE, "kz_tasks_check.cpp"), os.path.join(CSRC, "kz_tasks.hpp"),
            os.path.join(CSRC, "fft_core.hpp"), os.path.join(HERE, "hip", "hip_runtime.h")]
    if not os.path.exists(exe) or any(os.path.getmtime(s) > os.path.getmtime(exe) for s in srcs):
        cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
               "-I" + HERE, "-I" + CSRC, srcs[0], "-o", exe + ".tmp"]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, "compile failed:\n" + r.stdout[-3000:]
        os.replace(exe + ".tmp", exe)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout[-3000:]
