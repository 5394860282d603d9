"""Build the library's sources for the CPU emulation of HIP (tests only):
g++ with AddressSanitizer, the HIP shim of this folder in place of the HIP
headers.  Output: tests/cpuemu/_build/libgmg_emu.so."""
import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1904_03317_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libgmg_emu.so")
FLAGS = ["-std=c++20", "-O1", "-g", "-fPIC", "-pthread", "-fsanitize=address", "-fno-omit-frame-pointer",
         "-Wno-unknown-pragmas", "-Wno-unused-function", f"-I{HERE}", f"-I{ROOT}/include"]


def sources():
    host = [os.path.join(CSRC, "host", f) for f in sorted(os.listdir(os.path.join(CSRC, "host"))) if f.endswith(".cpp")]
    # mark.hip sorts with the device radix sort of hipcub; the emulation
    # takes mark_emu.cpp (same contract, a host sort) in its place
    dev = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip") and f != "mark.hip"]
    return host + dev + [os.path.join(HERE, "mark_emu.cpp")]


def _cc(src):
    obj = os.path.join(OUT, os.path.basename(os.path.dirname(src)) + "_" + os.path.basename(src) + ".o")
    cmd = ["g++", *FLAGS, "-x", "c++", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(" ".join(cmd) + "\n" + r.stderr[-4000:])
    return obj


def build(jobs=8):
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_cc, sources()))
    cmd = ["g++", "-shared", "-fsanitize=address", "-pthread", *objs, "-o", LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr[-4000:])
    return LIB


if __name__ == "__main__":
    print(build())
